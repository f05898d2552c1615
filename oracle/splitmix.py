"""SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) used as a counter-based generator.

The paper does not say how the ALS start tensor of a row absorption is
chosen; here it is filled with a deterministic pseudo-random tensor so that
the oracle and the GPU path start from the same point.  Both sides implement
the generator from its published definition:

    gamma = 0x9E3779B97F4A7C15
    mix(z): z = (z ^ z>>30) * 0xBF58476D1CE4E5B9
            z = (z ^ z>>27) * 0x94D049BB133111EB
            return z ^ z>>31
    n-th output of the stream with state s:  mix(s + (n+1)*gamma)   (mod 2^64)

A stream q of a run seeded with ``seed`` has state s_q = mix(seed + (q+1)*gamma);
its e-th value is mapped to [-1, 1) as  2*((x >> 11) * 2^-53) - 1.
"""
import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK = (1 << 64) - 1


def mix(z):
    """SplitMix64 output function on Python ints (exact mod 2^64)."""
    z &= MASK
    z = ((z ^ (z >> 30)) * M1) & MASK
    z = ((z ^ (z >> 27)) * M2) & MASK
    return z ^ (z >> 31)


def stream_state(seed, q):
    return mix(seed + (q + 1) * GAMMA)


def _mix_u64(z):
    # vectorised form of ``mix`` on uint64 arrays (wrapping arithmetic)
    z = z ^ (z >> np.uint64(30))
    z = z * np.uint64(M1)
    z = z ^ (z >> np.uint64(27))
    z = z * np.uint64(M2)
    return z ^ (z >> np.uint64(31))


def uniform(seed, q, count):
    """``count`` values in [-1, 1) from stream ``q``."""
    s = np.uint64(stream_state(seed, q))
    n = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = _mix_u64(s + n * np.uint64(GAMMA))
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0


def als_stream(side, row, col):
    """Stream id of the ALS start tensor for (side, absorbed row, column)."""
    return (side << 40) | (row << 20) | col
