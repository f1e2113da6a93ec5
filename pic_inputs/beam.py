"""Cold relativistic beam loader (the uniform drifting beam of Sec. 3).

Positions are stratified: every cell receives `ppc` points drawn uniformly
inside it, cells enumerated x-fastest, so particle p lives in cell p // ppc.
Momenta (u = gamma*v, per unit mass, c = 1) are u0 * (z_hat + sigma * xi)
with xi ~ N(0, I_3) and u0 = sqrt(gamma^2 - 1).  The beam axis is z.

Arrays are float64.  Layout: x has shape (N, dims) holding absolute positions
(2D: columns x, z; 3D: columns x, y, z), u has shape (N, 3) holding (ux, uy, uz).
"""
import numpy as np


def beam_weight(n0, cell_volume, ppc):
    """Macro-particle weight so that ppc particles per cell carry density n0."""
    return float(n0) * float(cell_volume) / float(ppc)


def load_beam(dims, n, ppc, gamma, sigma, seed, d=(1.0, 1.0, 1.0), cells=None):
    """Return (x, u) for a uniform beam on a periodic box.

    dims  : 2 or 3
    n     : (nx, nz) for 2D or (nx, ny, nz) for 3D cell counts
    ppc   : particles per cell
    gamma : beam Lorentz factor
    sigma : relative Gaussian momentum spread (applied to all 3 components)
    seed  : PCG64 seed
    d     : (dx, dz) or (dx, dy, dz) cell sizes
    cells : optional array of linear cell indices to load (default: all cells);
            lets a caller build a clumped or partial beam for edge cases.
    """
    n = tuple(int(v) for v in n)
    d = tuple(float(v) for v in d)
    assert dims in (2, 3) and len(n) == dims and len(d) >= dims
    rng = np.random.Generator(np.random.PCG64(seed))
    ncell = int(np.prod(n))
    if cells is None:
        cells = np.arange(ncell, dtype=np.int64)
    cells = np.asarray(cells, dtype=np.int64)
    npart = cells.size * ppc
    cid = np.repeat(cells, ppc)
    # decompose linear cell index, x fastest
    coords = []
    rem = cid
    for a in range(dims):
        coords.append(rem % n[a])
        rem = rem // n[a]
    r = rng.random((npart, dims))
    x = np.empty((npart, dims), dtype=np.float64)
    for a in range(dims):
        x[:, a] = (coords[a] + r[:, a]) * d[a]
    u0 = np.sqrt(gamma * gamma - 1.0)
    xi = rng.standard_normal((npart, 3))
    u = np.empty((npart, 3), dtype=np.float64)
    u[:, 0] = u0 * sigma * xi[:, 0]
    u[:, 1] = u0 * sigma * xi[:, 1]
    u[:, 2] = u0 * (1.0 + sigma * xi[:, 2])
    return x, u
