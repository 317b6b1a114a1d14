"""The oracle on small periodic windows of a large lattice.

One time step changes a site's distributions through its neighbours' lapse
and metric (the derivative stencil) and through streaming, so information
moves at most two sites per step (Chebyshev distance), and the output moments
reach one site further (their half-source uses the stencil once more); the
initialisation from fields uses the stencil once.  So after `steps` steps from
fields, the moments and distributions at the centre of a periodic window of
radius R = 2 * steps + 2 cut from the initial fields are those of the whole
lattice at that site: the window's own wrap-around reaches the centre only
later.  This gives exact oracle values at sampled sites of lattices far too
large for the oracle to evolve whole.
"""

import numpy as np

import oracle


def window_radius(steps: int) -> int:
    return 2 * steps + 2


def cut(u: np.ndarray, centre, R: int) -> np.ndarray:
    """The fields u[:, z-R..z+R, y-R..y+R, x-R..x+R] with periodic wrap."""
    nz, ny, nx = u.shape[1:]
    z, y, x = centre
    iz = np.arange(z - R, z + R + 1) % nz
    iy = np.arange(y - R, y + R + 1) % ny
    ix = np.arange(x - R, x + R + 1) % nx
    return np.ascontiguousarray(u[np.ix_(np.arange(u.shape[0]), iz, iy, ix)])


def sampled(u0: np.ndarray, centres, tau: float, steps: int, slicing=oracle.HARMONIC,
            collision=oracle.COLLISION_BGK, R: int | None = None):
    """Oracle moments (16, S) and distributions (16, 19, S) at `centres`
    ((z, y, x) triples) after `steps` steps of the D3Q19 step from u0."""
    R = window_radius(steps) if R is None else R
    w = 2 * R + 1
    us, fs = [], []
    for c in centres:
        o = oracle.Oracle(w, w, w, tau, slicing, collision=collision)
        o.init_fields(cut(u0, c, R))
        o.step(steps)
        us.append(o.moments()[:, R, R, R])
        fs.append(o.distributions()[:, :, R, R, R])
        o.close()
    return np.stack(us, axis=-1), np.stack(fs, axis=-1)


def sample_centres(n: int, count: int, seed: int):
    """Corner and face sites of an n^3 lattice (where the periodic wrap acts)
    and `count` seeded random sites, as (z, y, x) triples."""
    rng = np.random.Generator(np.random.PCG64(seed))
    edge = [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, n // 2), (n - 1, 0, 1), (n // 2, n // 2, 0),
            (1, n - 2, n - 1)]
    return edge + [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(count)]
