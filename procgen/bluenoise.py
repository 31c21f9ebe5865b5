"""Blue-noise threshold texture by void-and-cluster (Ulichney, "The void-and-cluster method for
dither array generation", SPIE 1993), written from the published description.

The texture is a table of the random numbers the sampling step draws (one threshold per
pixel, tiled over the frame), so it is an input like the scene: both the GPU path and the
oracle take it as given.  Energies are integer sums of a quantised toroidal Gaussian, so the
result does not depend on summation order; ties go to the lowest linear index.
"""
import numpy as np


def _kernel(T: int, sigma: float):
    d = np.minimum(np.arange(T), T - np.arange(T)).astype(np.float64)
    g = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2.0 * sigma * sigma))
    return np.round(g * (1 << 20)).astype(np.int64)


def void_and_cluster(T: int = 64, sigma: float = 1.5, seed: int = 0, init_frac: float = 0.1):
    """Rank matrix [T, T] (a permutation of 0 .. T*T-1): thresholding at rank < m gives a
    well-spread pattern of m pixels for every m."""
    K = _kernel(T, sigma)
    flatK = K.reshape(-1)

    def splat(E, i, sgn):
        y, x = divmod(int(i), T)
        E += sgn * np.roll(np.roll(K, y, 0), x, 1)

    rng = np.random.default_rng([int(seed), 0xB1E])
    n1 = max(1, int(init_frac * T * T))
    B = np.zeros((T, T), bool)
    B.flat[rng.choice(T * T, n1, replace=False)] = True
    E = np.zeros((T, T), np.int64)
    for i in np.flatnonzero(B):
        splat(E, i, 1)
    lo, hi = np.iinfo(np.int64).min, np.iinfo(np.int64).max
    tightest = lambda B, E: int(np.argmax(np.where(B, E, lo)))     # 1 with the most 1-energy
    largest_void = lambda B, E: int(np.argmin(np.where(B, hi, E)))  # 0 with the least 1-energy
    # initial pattern: move the tightest cluster into the largest void until they coincide
    for _ in range(T * T):
        c = tightest(B, E)
        B.flat[c] = False
        splat(E, c, -1)
        v = largest_void(B, E)
        B.flat[v] = True
        splat(E, v, 1)
        if v == c:
            break
    rank = np.full(T * T, -1, np.int64)
    # phase 1: remove the initial points tightest-first, ranks n1-1 .. 0
    B1, E1 = B.copy(), E.copy()
    for r in range(n1 - 1, -1, -1):
        c = tightest(B1, E1)
        rank[c] = r
        B1.flat[c] = False
        splat(E1, c, -1)
    # phases 2 and 3: fill the largest void, ranks n1 .. T*T-1 (with a linear energy the
    # tightest cluster of 0s is the 0 with the least 1-energy, so phase 3 is the same rule)
    B2, E2 = B.copy(), E.copy()
    for r in range(n1, T * T):
        v = largest_void(B2, E2)
        rank[v] = r
        B2.flat[v] = True
        splat(E2, v, 1)
    assert (rank >= 0).all()
    return rank.reshape(T, T)


def blue_noise_thresholds(T: int = 64, seed: int = 0):
    """float32 [T, T] thresholds u = (rank + 1/2) / T^2 in (0, 1), exact in binary32."""
    return ((void_and_cluster(T, seed=seed).astype(np.float64) + 0.5) / (T * T)).astype(np.float32)
