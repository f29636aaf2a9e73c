"""SplitMix64 as a counter-based generator (oracle side).

Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014: a generator with seed ``s`` returns ``mix64(s + k * GAMMA)`` for
k = 1, 2, ...; ``mix64`` is their variant-13 finaliser.  Output ``n`` (0-based)
of the stream with seed ``s`` is therefore ``mix64(s + (n + 1) * GAMMA)``.

Ray jitter: for box key b, cast axis w, cell (i, j) the counter is
``n = 2 * ((b << 32) | (w << 30) | (i << 15) | j) + c`` with c = 0 for the u
jitter and c = 1 for the v jitter; the jitter is the top 24 bits times 2^-24
(exact in float32 and float64).
"""
import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK = (1 << 64) - 1


def mix64(z):
    """Variant-13 finaliser on Python ints (reference scalar form)."""
    z &= MASK
    z = ((z ^ (z >> 30)) * M1) & MASK
    z = ((z ^ (z >> 27)) * M2) & MASK
    return z ^ (z >> 31)


def splitmix64(seed, n):
    """Output n (0-based) of the SplitMix64 stream with the given seed (scalar)."""
    return mix64((seed + (n + 1) * GAMMA) & MASK)


def splitmix64_np(seed, n):
    """Vectorised splitmix64 over a uint64 array of counters (wrap-around arithmetic)."""
    n = np.asarray(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK) + (n + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        z = z ^ (z >> np.uint64(31))
    return z


def u24(x):
    """Top 24 bits of a uint64 as a float64 in [0, 1)."""
    return (np.asarray(x, dtype=np.uint64) >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)


def ray_counter(box_key, w, i, j):
    i = np.asarray(i, dtype=np.uint64)
    j = np.asarray(j, dtype=np.uint64)
    return ((np.uint64(box_key) << np.uint64(32)) | (np.uint64(w) << np.uint64(30))
            | (i << np.uint64(15)) | j)


def jitter(seed, box_key, w, i, j):
    """(xi, eta) in [0,1)^2 for the cells (i, j) of cast axis w of box ``box_key``."""
    key = ray_counter(box_key, w, i, j)
    with np.errstate(over="ignore"):
        xi = u24(splitmix64_np(seed, np.uint64(2) * key))
        eta = u24(splitmix64_np(seed, np.uint64(2) * key + np.uint64(1)))
    return xi, eta
