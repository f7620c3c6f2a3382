"""Counter-based SplitMix64 (Steele, Lea and Flood, 2014) for seeded inputs.

Output k of the stream seeded with s is mix(s + (k + 1) * 0x9E3779B97F4A7C15)
with mix the SplitMix64 finaliser; the uniform variate on [-1, 1) takes the
top 53 bits.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, counter):
    """Vectorised k-th output (k = counter) of the stream seeded with seed."""
    with np.errstate(over="ignore"):
        k = np.asarray(counter, dtype=np.uint64)
        z = np.uint64(seed) + (k + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        return z ^ (z >> np.uint64(31))


def uniform_pm1(seed, counter):
    z = splitmix64(seed, counter)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0


def perturbation(shape, seed, amplitude, solid=None):
    """Velocity field [3][nz][ny][nx]: amplitude * xi, xi ~ U[-1,1) from
    counter 3*cell + component; zero in solid cells."""
    nx, ny, nz = shape
    N = nx * ny * nz
    cell = np.arange(N, dtype=np.uint64)
    u = np.empty((3, N))
    for d in range(3):
        u[d] = amplitude * uniform_pm1(seed, np.uint64(3) * cell + np.uint64(d))
    if solid is not None:
        u[:, np.asarray(solid).reshape(-1).astype(bool)] = 0.0
    return u.reshape(3, nz, ny, nx)
