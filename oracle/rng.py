"""Counter-based normal draws used by the method (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method draws random numbers in two places: the Gaussian test matrix of the
HMT range finder in the initialisation, and the random perturbation xi_t of the
rank safeguard (supplement, "Initialization" and "Ensuring Sufficient Precision
in the Proximal Operation").  Both sides of the parity test implement the same
published generator independently, so the draws agree:

* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): state x advances by the golden
  gamma 0x9E3779B97F4A7C15 and each output is the state passed through the
  variant-13 finaliser mix64.
* For a (seed, stream) pair the start state is
  x0 = seed XOR (stream * 0xD1B54A32D192ED03)  (mod 2^64);
  draw number c (c = 0, 1, ...) is mix64(x0 + (c + 1) * gamma).
* A uniform in (0, 1) is ((v >> 11) + 0.5) * 2^-53.
* Normal number i is Box-Muller on draws 2i and 2i+1:
  sqrt(-2 ln u1) * cos(2 pi u2).
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_SKEW = np.uint64(0xD1B54A32D192ED03)

STREAM_SKETCH = 1          # HMT test matrix, entry (i, j) of an m x k0 matrix -> index i*k0 + j
STREAM_SAFEGUARD = 0x100   # + outer iteration t; entry i of an m-vector -> index i


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def raw_draws(seed: int, stream: int, count: int) -> np.ndarray:
    """The 64-bit outputs: draw c is mix64(x0 + (c + 1) * gamma)."""
    with np.errstate(over="ignore"):
        x0 = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ (np.uint64(stream & 0xFFFFFFFFFFFFFFFF) * _SKEW)
        c = np.arange(1, count + 1, dtype=np.uint64)
        return _mix64(x0 + c * _GAMMA)


def uniform_draws(seed: int, stream: int, count: int) -> np.ndarray:
    v = raw_draws(seed, stream, count)
    return ((v >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def normals(seed: int, stream: int, count: int) -> np.ndarray:
    u = uniform_draws(seed, stream, 2 * count)
    u1, u2 = u[0::2], u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
