"""Counter-based SplitMix64 stream (Steele, Lea and Flood, OOPSLA 2014).

Every random draw used to build a workload comes from here, so a seed fully
determines a mesh and its initial data on any machine.
"""

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, start: int, n: int) -> np.ndarray:
    """Outputs number start..start+n-1 of the SplitMix64 sequence seeded by `seed`."""
    with np.errstate(over="ignore"):
        ctr = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + ctr * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


class Stream:
    """Sequential view of one SplitMix64 sequence."""

    def __init__(self, seed: int):
        self.seed = int(seed)
        self.pos = 0

    def bits(self, n: int) -> np.ndarray:
        out = splitmix64(self.seed, self.pos, n)
        self.pos += n
        return out

    def uniform(self, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        """n doubles uniform in [lo, hi): top 53 bits scaled by 2^-53."""
        u = (self.bits(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        return lo + (hi - lo) * u

    def log_uniform(self, n: int, lo: float, hi: float) -> np.ndarray:
        return np.exp(self.uniform(n, np.log(lo), np.log(hi)))
