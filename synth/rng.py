"""Counter-based SplitMix64 streams (Steele, Lea & Flood 2014; the mixing
constants are those of the published SplitMix64 finaliser).

Value k (k = 0, 1, ...) of the stream with seed ``s`` is the (k+1)-th output
of a sequential SplitMix64 started from state ``s``, so a stream can be drawn
in any order or in bulk.  Uniforms use the top 53 bits; normals use
Box-Muller on pairs of uniforms.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

BASE_SEED = 1805021440


def _mix(z):
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_seed(seed, stream_id):
    """Sub-stream seed = seed xor (stream_id * GAMMA) (mod 2**64)."""
    with np.errstate(over="ignore"):
        return np.uint64(seed) ^ (np.uint64(stream_id) * GAMMA)


class Stream:
    def __init__(self, seed, stream_id=0):
        self.state = stream_seed(seed, stream_id)
        self.k = 0

    def u64(self, n):
        with np.errstate(over="ignore"):
            idx = np.arange(self.k + 1, self.k + 1 + n, dtype=np.uint64)
            out = _mix(self.state + idx * GAMMA)
        self.k += n
        return out

    def uniform(self, n):
        return (self.u64(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def normal(self, n):
        m = (n + 1) // 2
        u1 = self.uniform(m)
        u2 = self.uniform(m)
        u1 = np.where(u1 <= 0.0, 2.0 ** -53, u1)
        r = np.sqrt(-2.0 * np.log(u1))
        z = np.concatenate([r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)])
        return z[:n]

    def integers(self, n, high):
        """Uniform integers in [0, high) (multiply-shift on 53-bit uniforms)."""
        return np.floor(self.uniform(n) * high).astype(np.int64)
