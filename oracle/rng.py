"""SplitMix64 counter-based generator — oracle side (test infrastructure only).

The method draws random sample positions (Alg. 2, first step: "pick a random
set of samples").  To make the GPU library and the oracle draw the SAME
positions without sharing code, each side implements the published SplitMix64
generator (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; the constants are those of S. Vigna's public
``splitmix64.c``) in counter form:

    value(seed, c) = mix(seed + (c + 1) * GAMMA)   (mod 2**64)

which is the (c+1)-th output of a SplitMix64 stream started from state ``seed``.

Counter layout (a reading of the paper, which does not fix the distribution):

* random samples of bond b in sweep s, sample j:  c = s * 2**40 + b * 2**24 + j
* rank-1 start, sample q, mode k:                 c = 2**63 + q * 2**16 + k
* Monte Carlo estimator j, point i, coordinate k (m coordinates per point):
                                                  c = 2**62 + j * 2**40 + i * m + k
* lattice shift of estimator j, coordinate k:     c = 2**62 + 2**61 + j * 2**6 + k

A uniform integer in [0, N), N < 2**32, is ``((u >> 32) * N) >> 32``; a
uniform double in the open interval (0, 1) is ``((u >> 11) + 0.5) * 2**-53``.

Pinned by: the published first outputs of the seed-0 stream (tests/golden).
"""

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB

START_DOMAIN = 1 << 63


def mix(z):
    """SplitMix64 output function applied to a 64-bit state."""
    z &= MASK
    z = ((z ^ (z >> 30)) * M1) & MASK
    z = ((z ^ (z >> 27)) * M2) & MASK
    return z ^ (z >> 31)


def value(seed, counter):
    """(counter+1)-th output of the SplitMix64 stream whose state starts at seed."""
    return mix((seed + ((counter + 1) * GAMMA)) & MASK)


def stream(seed, count):
    """First ``count`` outputs of the sequential SplitMix64 stream (for pins)."""
    x = seed & MASK
    out = []
    for _ in range(count):
        x = (x + GAMMA) & MASK
        out.append(mix(x))
    return out


def uniform_index(u, n):
    """Map a 64-bit draw to [0, n) with the high 32 bits (n < 2**32)."""
    assert 0 < n < (1 << 32)
    return ((u >> 32) * n) >> 32


def sample_counter(sweep, bond, j):
    return (sweep << 40) + (bond << 24) + j


def start_counter(q, k):
    return START_DOMAIN + (q << 16) + k


MC_DOMAIN = 1 << 62
SHIFT_DOMAIN = (1 << 62) + (1 << 61)


def mc_counter(j, i, m, k):
    return MC_DOMAIN + (j << 40) + i * m + k


def shift_counter(j, k):
    return SHIFT_DOMAIN + (j << 6) + k


def uniform_open01(u):
    """A 64-bit draw mapped to a double in (0, 1): the top 53 bits, centred in their cell."""
    return ((u >> 11) + 0.5) * 2.0 ** -53
