"""SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) -- the oracle's own implementation.

The solver draws one vector q_j per greedy step j to build its initial ALS
vector (the paper leaves the choice open in Algorithm 1: "pick initial
vector v").  Stream ``j`` of seed ``s`` starts from the state
s XOR (j * 0xD1B54A32D192ED03) mod 2^64; output k >= 1 is the SplitMix64
finaliser applied to state + k * 0x9E3779B97F4A7C15, and its top 53 bits
map to a double in [-1, 1) as (z >> 11) * 2^-52 - 1.
"""
import numpy as np

GOLDEN_GAMMA = 0x9E3779B97F4A7C15
STREAM_MUL = 0xD1B54A32D192ED03
_M64 = (1 << 64) - 1


def mix64(z: int) -> int:
    """The SplitMix64 output finaliser on a Python int (mod 2^64)."""
    z &= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def splitmix64_sequence(state: int, n: int):
    """First n outputs of SplitMix64 started from ``state`` (Python ints)."""
    out = []
    for k in range(1, n + 1):
        out.append(mix64(state + k * GOLDEN_GAMMA))
    return out


def uniform_pm1(seed: int, stream: int, n: int) -> np.ndarray:
    """n doubles in [-1, 1) from stream ``stream`` of ``seed`` (vectorised)."""
    state = (int(seed) ^ ((int(stream) * STREAM_MUL) & _M64)) & _M64
    k = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(state) + k * np.uint64(GOLDEN_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0
