"""Counter-based splitmix64 streams in numpy uint64 arithmetic.

splitmix64 (Steele, Lea, Flood, OOPSLA 2014): state advances by the golden
gamma 0x9E3779B97F4A7C15 and each output is the state passed through the
variant-13 finaliser (shifts 30/27/31, multipliers 0xBF58476D1CE4E5B9 and
0x94D049BB133111EB).  Element i of a stream is the finaliser applied to
base + (i + 1) * gamma, so any slice of a stream can be produced directly.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    """The splitmix64 finaliser, elementwise on a uint64 array (wrapping)."""
    z = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def _base(seed, stream):
    with np.errstate(over="ignore"):
        s = splitmix64(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))
        t = splitmix64(np.array([(stream * 0x632BE59BD9B4E019) & 0xFFFFFFFFFFFFFFFF],
                                dtype=np.uint64))
        return splitmix64(s ^ t)[0]


def stream_u64(seed, stream, count, start=0):
    """Elements [start, start+count) of the splitmix64 stream (seed, stream)."""
    base = _base(seed, stream)
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return splitmix64(base + idx * _GAMMA)


def stream_uniform(seed, stream, count, start=0):
    """Uniform doubles in [0, 1) from the top 53 bits of the u64 stream."""
    u = stream_u64(seed, stream, count, start)
    return (u >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
